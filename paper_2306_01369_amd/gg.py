"""Thin Python binding of libgg (include/gg.h): argument marshalling only.

Every step of the simulation runs in the HIP kernels behind the C ABI; this
module converts NumPy arrays / torch tensors to pointers and status codes to
exceptions.  It fails loudly when the library has not been built: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgg.so")

GG_OK, GG_ERR_INVALID, GG_ERR_OOM, GG_ERR_HIP, GG_ERR_CAPACITY, GG_ERR_NONFINITE, GG_ERR_NO_TAPE, \
    GG_ERR_UNSUPPORTED = range(8)
GG_MEM_HOST, GG_MEM_DEVICE = 0, 1
GG_FLAG_PROFILE, GG_FLAG_DIAGNOSTICS, GG_FLAG_TAPE, GG_FLAG_GRAPH, GG_FLAG_FUSED = 1, 2, 4, 8, 16
FIELD = {"pos": 0, "vel": 1, "cell_index": 2, "contacts": 3, "impulses": 4, "stats": 5, "dv": 6,
         "radius": 7, "body_poses": 8}
SHAPES = {"plane": 0, "box": 1, "capsule": 2, "grid": 3}

EXPORTS = ("gg_create", "gg_set_bodies", "gg_set_grids", "gg_step", "gg_step_backward", "gg_read",
           "gg_render_depth", "gg_goal_reward", "gg_goal_reward_noalloc", "gg_destroy",
           "gg_status_string", "gg_error_detail")


class GGError(RuntimeError):
    def __init__(self, status, detail):
        self.status = status
        super().__init__(f"gg status {status}: {detail}")


class CapacityError(GGError):
    pass


class Body(C.Structure):
    _fields_ = [("env", C.c_int32), ("shape", C.c_int32), ("params", C.c_float * 4),
                ("pose", C.c_float * 12), ("twist", C.c_float * 6)]


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("origin", C.c_float * 3),
                ("inv_spacing", C.c_float), ("offset", C.c_int64)]


class Camera(C.Structure):
    _fields_ = [("env", C.c_int32), ("kind", C.c_int32), ("width", C.c_int32), ("height", C.c_int32),
                ("pose", C.c_float * 12), ("params", C.c_float * 4)]


CAMERA_KINDS = {"ortho": 0, "perspective": 1}


def make_cameras(cams):
    """gg_camera array from dicts {"env", "kind" ("ortho" | "perspective"),
    "width", "height", "pose" (3 x 4, camera -> world), "params" (p0, p1, far)}."""
    arr = (Camera * max(1, len(cams)))()
    for k, c in enumerate(cams):
        A = arr[k]
        A.env = int(c.get("env", 0))
        A.kind = CAMERA_KINDS[c["kind"]] if isinstance(c["kind"], str) else int(c["kind"])
        A.width, A.height = int(c["width"]), int(c["height"])
        pose = np.asarray(c["pose"], np.float64).reshape(12)
        for q in range(12):
            A.pose[q] = float(pose[q])
        prm = list(c["params"]) + [0.0] * (4 - len(c["params"]))
        for q in range(4):
            A.params[q] = float(prm[q])
    return arr


class Params(C.Structure):
    _fields_ = [("dt", C.c_float), ("alpha", C.c_float), ("mu", C.c_float), ("gravity", C.c_float * 3),
                ("n_iters", C.c_int32), ("cell_size", C.c_float), ("hash_size", C.c_int64),
                ("relax", C.c_float), ("mass_split", C.c_int32), ("checkpoint_every", C.c_int32),
                ("max_contacts_per_particle", C.c_int32), ("precision", C.c_int32),
                ("density", C.c_float), ("flags", C.c_uint32), ("reorder_every", C.c_int32),
                ("tile_max_cells", C.c_int32), ("tile_max_stage", C.c_int32),
                ("tile_node_shift", C.c_int32), ("tile_threads", C.c_int32), ("cyclic_z", C.c_float * 2),
                ("pja_lanes", C.c_int32), ("device", C.c_int32),
                ("stream", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("steps_done", C.c_int64), ("steps_total", C.c_int64), ("n_pp", C.c_int64),
                ("n_pb", C.c_int64), ("candidates", C.c_int64), ("max_contacts", C.c_int64),
                ("capacity", C.c_int64), ("last_status", C.c_int64), ("n", C.c_int64),
                ("n_buckets", C.c_int64), ("ms_detect", C.c_double), ("ms_pja", C.c_double),
                ("ms_integrate", C.c_double), ("pja_launches", C.c_int64),
                ("contacts_summed", C.c_int64), ("detect_fallback", C.c_int64),
                ("detect_items", C.c_int64), ("device_bytes_peak", C.c_int64),
                ("tile_threads", C.c_int32), ("tile_node_shift", C.c_int32), ("tile_max_cells", C.c_int32),
                ("tile_max_stage", C.c_int32), ("detect_workgroups", C.c_int32), ("reorder_every", C.c_int32),
                ("pja_lanes", C.c_int32), ("detect_queues", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_LIB = None


def lib():
    """Load libgg.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(there is no CPU fallback)")
        # torch bundles its own HIP runtime with the same soname; load it first so
        # that a process using both shares one runtime (two runtimes in one
        # process cannot both open the device).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.gg_create.restype = i32
        L.gg_create.argtypes = [C.POINTER(Params), i32, vp, i64, vp, vp, vp, i32, C.POINTER(vp)]
        L.gg_set_bodies.restype = i32
        L.gg_set_bodies.argtypes = [vp, i32, vp, i32]
        L.gg_set_grids.restype = i32
        L.gg_set_grids.argtypes = [vp, i32, vp, i64, vp, i32]
        L.gg_step.restype = i32
        L.gg_step.argtypes = [vp, i32, vp, i32]
        L.gg_step_backward.restype = i32
        L.gg_step_backward.argtypes = [vp, vp, vp, vp, vp, vp, i32]
        L.gg_read.restype = i32
        L.gg_read.argtypes = [vp, i32, vp, i64, C.POINTER(i64), i32]
        L.gg_render_depth.restype = i32
        L.gg_render_depth.argtypes = [vp, i32, vp, vp, i64, i32]
        L.gg_goal_reward.restype = i32
        L.gg_goal_reward.argtypes = [vp, vp, vp, vp, i32]
        L.gg_goal_reward_noalloc.restype = i32
        L.gg_goal_reward_noalloc.argtypes = [vp, vp, vp, vp, i32]
        L.gg_destroy.restype = None
        L.gg_destroy.argtypes = [vp]
        L.gg_status_string.restype = C.c_char_p
        L.gg_status_string.argtypes = [i32]
        L.gg_error_detail.restype = C.c_char_p
        L.gg_error_detail.argtypes = []
        _LIB = L
    return _LIB


def _check(st):
    if st != GG_OK:
        detail = lib().gg_error_detail().decode()
        if st == GG_ERR_CAPACITY:
            raise CapacityError(st, detail)
        raise GGError(st, detail)


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _arg(a, dtype, shape=None):
    """(pointer, where, keepalive) for a NumPy array or a torch tensor."""
    if a is None:
        return None, GG_MEM_HOST, None
    if _is_torch(a):
        import torch
        tdt = {np.float32: torch.float32, np.int64: torch.int64}[dtype]
        t = a.detach()
        if t.dtype != tdt:
            t = t.to(tdt)
        t = t.contiguous()
        return C.c_void_p(t.data_ptr()), (GG_MEM_DEVICE if t.is_cuda else GG_MEM_HOST), t
    arr = np.ascontiguousarray(np.asarray(a, dtype=dtype))
    if shape is not None:
        arr = arr.reshape(shape)
    return arr.ctypes.data_as(C.c_void_p), GG_MEM_HOST, arr


def make_body(d):
    """gg_body from a scenes-style dict (shape, params, R, t, nu, omega, env)."""
    b = Body()
    b.env = int(d.get("env", 0))
    b.shape = SHAPES[d["shape"]] if isinstance(d["shape"], str) else int(d["shape"])
    for q in range(4):
        b.params[q] = float(d["params"][q])
    R = np.asarray(d["R"], np.float64).reshape(3, 3)
    t = np.asarray(d["t"], np.float64)
    for r in range(3):
        for c in range(3):
            b.pose[4 * r + c] = float(R[r, c])
        b.pose[4 * r + 3] = float(t[r])
    for q in range(3):
        b.twist[q] = float(d["nu"][q])
        b.twist[3 + q] = float(d["omega"][q])
    return b


class Sim:
    """One gg_sim handle.  Positions/velocities/radii may be NumPy arrays (host)
    or torch tensors (host or device)."""

    def __init__(self, x, v, radius, bodies=(), *, dt=1e-3, alpha=0.2, mu=0.5, n_iters=20,
                 gravity=(0.0, 0.0, -9.81), cell_size=0.0, hash_size=0, relax=1.0, mass_split=True,
                 max_contacts=0, density=2500.0, env_offsets=None, device=0, stream=None,
                 profile=False, diagnostics=False, reorder_every=0, tile_max_cells=0,
                 tile_max_stage=0, tile_node_shift=0, tile_threads=0, differentiable=False, checkpoint_every=0,
                 graph=False, precision=0, cyclic_z=None, fused=False, pja_lanes=0):
        L = lib()
        P = Params()
        P.dt, P.alpha, P.mu = dt, alpha, mu
        for a in range(3):
            P.gravity[a] = gravity[a]
        P.n_iters = n_iters
        P.cell_size = cell_size
        P.hash_size = int(hash_size)
        P.relax = relax
        P.mass_split = 1 if mass_split else 0
        P.max_contacts_per_particle = int(max_contacts)
        P.density = density
        P.flags = (GG_FLAG_PROFILE if profile else 0) | (GG_FLAG_DIAGNOSTICS if diagnostics else 0) | \
            (GG_FLAG_TAPE if differentiable else 0) | (GG_FLAG_GRAPH if graph else 0) | \
            (GG_FLAG_FUSED if fused else 0)
        P.checkpoint_every = int(checkpoint_every)
        P.precision = int(precision)
        P.reorder_every = int(reorder_every)
        P.tile_max_cells = int(tile_max_cells)
        P.tile_max_stage = int(tile_max_stage)
        P.tile_node_shift = int(tile_node_shift)
        P.tile_threads = int(tile_threads)
        P.pja_lanes = int(pja_lanes)
        if cyclic_z is not None:
            P.cyclic_z[0], P.cyclic_z[1] = float(cyclic_z[0]), float(cyclic_z[1])
        P.device = device
        P.stream = stream
        n = int(x.shape[0])
        px, wx, kx = _arg(x, np.float32, (-1, 3))
        pv, wv, kv = _arg(v, np.float32, (-1, 3))
        pr, wr, kr = _arg(radius, np.float32)
        if len({wx, wv, wr}) != 1:
            raise ValueError("x, v and radius must all live on the host or all on the device")
        offs = None
        n_envs = 1
        if env_offsets is not None:
            offs = np.ascontiguousarray(env_offsets, np.int64)
            n_envs = len(offs) - 1
        h = C.c_void_p()
        st = L.gg_create(C.byref(P), n_envs, None if offs is None else offs.ctypes.data_as(C.c_void_p), n,
                         px, pv, pr, wx, C.byref(h))
        _check(st)
        self._h = h
        self.n = n
        self.n_envs = n_envs
        self.params = P
        self.n_bodies = 0
        if bodies:
            self.set_bodies(bodies)

    def close(self):
        if getattr(self, "_h", None):
            lib().gg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_bodies(self, bodies):
        """Bodies as scenes-style dicts (or gg_body records).  A "grid" body
        carries its samples: d["grid"] = {"values": (nz, ny, nx) float32,
        "origin": (3,), "inv_spacing": float}; the distinct grids are
        registered (gg_set_grids) and indexed through params[0]."""
        bodies = list(bodies)
        grids, index, recs = [], {}, []
        for b in bodies:
            if isinstance(b, dict) and b.get("shape") == "grid":
                g = b["grid"]
                key = id(g["values"])
                if key not in index:
                    index[key] = len(grids)
                    grids.append(g)
                b = dict(b, params=[float(index[key]), 0.0, 0.0, 0.0])
            recs.append(make_body(b) if isinstance(b, dict) else b)
        if grids:
            self.set_grids(grids)
        arr = (Body * max(1, len(recs)))(*recs)
        _check(lib().gg_set_bodies(self._h, len(recs), arr, GG_MEM_HOST))
        self.n_bodies = len(recs)

    def set_grids(self, grids):
        """Register SDF grids: list of {"values": (nz, ny, nx), "origin", "inv_spacing"}."""
        descs = (Grid * max(1, len(grids)))()
        chunks, off = [], 0
        for k, g in enumerate(grids):
            vals = np.ascontiguousarray(g["values"], np.float32)
            nz, ny, nx = vals.shape
            d = descs[k]
            d.nx, d.ny, d.nz = nx, ny, nz
            for a in range(3):
                d.origin[a] = float(g["origin"][a])
            d.inv_spacing = float(g["inv_spacing"])
            d.offset = off
            chunks.append(vals.ravel())
            off += vals.size
        allv = np.concatenate(chunks) if chunks else np.zeros(1, np.float32)
        _check(lib().gg_set_grids(self._h, len(grids), descs, int(off), allv.ctypes.data_as(C.c_void_p),
                                  GG_MEM_HOST))
        self._grids = list(grids)

    def step(self, n_steps=1, twists=None):
        if twists is not None:
            size = int(twists.numel()) if _is_torch(twists) else int(np.asarray(twists).size)
            if size != int(n_steps) * self.n_bodies * 6:
                raise ValueError(f"twists must hold n_steps x n_bodies x 6 = {int(n_steps)} x {self.n_bodies} x 6 "
                                 f"values, got {size}")
        pt, wt, kt = _arg(twists, np.float32)
        self.last_steps = int(n_steps)
        _check(lib().gg_step(self._h, int(n_steps), pt, wt))

    def read_bytes(self, field):
        w = C.c_int64(0)
        _check(lib().gg_read(self._h, FIELD[field], None, 0, C.byref(w), GG_MEM_HOST))
        return int(w.value)

    def read(self, field, out=None):
        """NumPy copy of a field, or copy into a given device tensor ``out``."""
        nbytes = self.read_bytes(field)
        if out is not None:
            w = C.c_int64(0)
            _check(lib().gg_read(self._h, FIELD[field], C.c_void_p(out.data_ptr()),
                                 out.numel() * out.element_size(), C.byref(w),
                                 GG_MEM_DEVICE if out.is_cuda else GG_MEM_HOST))
            return out
        if field == "stats":
            s = Stats()
            w = C.c_int64(0)
            _check(lib().gg_read(self._h, FIELD[field], C.byref(s), C.sizeof(s), C.byref(w), GG_MEM_HOST))
            return s.as_dict()
        dtype, cols = {"pos": (np.float32, 3), "vel": (np.float32, 3), "dv": (np.float32, 3),
                       "radius": (np.float32, 0), "cell_index": (np.int64, 0), "contacts": (np.int32, 2),
                       "impulses": (np.float32, 3), "body_poses": (np.float32, 12)}[field]
        item = np.dtype(dtype).itemsize * max(cols, 1)
        rows = nbytes // item
        arr = np.empty((rows, cols) if cols else (rows,), dtype)
        w = C.c_int64(0)
        if nbytes:
            _check(lib().gg_read(self._h, FIELD[field], arr.ctypes.data_as(C.c_void_p), nbytes, C.byref(w),
                                 GG_MEM_HOST))
        if field == "body_poses":
            return arr.reshape(-1, 3, 4)
        return arr

    def stats(self):
        return self.read("stats")

    def render_depth(self, cams, out=None):
        """Depth images of the current state (Sec. III-A observations): a list of
        (height, width) float32 arrays, or, with ``out`` (a device tensor of at
        least the total pixel count), the concatenated images written there."""
        A = make_cameras(cams)
        sizes = [int(c["width"]) * int(c["height"]) for c in cams]
        total = sum(sizes)
        if out is not None:
            _check(lib().gg_render_depth(self._h, len(cams), C.byref(A), C.c_void_p(out.data_ptr()),
                                         out.numel() * out.element_size(),
                                         GG_MEM_DEVICE if out.is_cuda else GG_MEM_HOST))
            return out
        buf = np.empty(total, np.float32)
        _check(lib().gg_render_depth(self._h, len(cams), C.byref(A), buf.ctypes.data_as(C.c_void_p), total * 4,
                                     GG_MEM_HOST))
        imgs, at = [], 0
        for c, m in zip(cams, sizes):
            imgs.append(buf[at:at + m].reshape(int(c["height"]), int(c["width"])))
            at += m
        return imgs

    def render_cameras(self, cam_array, n_cams, out):
        """Render a prepared gg_camera array (``make_cameras``) into ``out``, a
        float32 NumPy array or torch tensor (host or device) holding at least
        the total pixel count."""
        if _is_torch(out):
            ptr, nbytes = C.c_void_p(out.data_ptr()), out.numel() * out.element_size()
            where = GG_MEM_DEVICE if out.is_cuda else GG_MEM_HOST
        else:
            assert out.dtype == np.float32 and out.flags.c_contiguous
            ptr, nbytes, where = out.ctypes.data_as(C.c_void_p), out.nbytes, GG_MEM_HOST
        _check(lib().gg_render_depth(self._h, int(n_cams), C.byref(cam_array), ptr, nbytes, where))
        return out

    def goal_reward(self, boxes, noalloc=False):
        """(reward, inside) per environment for goal boxes n_envs x (lo, hi);
        noalloc: through gg_goal_reward_noalloc (no device allocation)."""
        bx = np.ascontiguousarray(boxes, np.float32).reshape(-1, 6)
        ne = bx.shape[0]
        if ne != self.n_envs:
            raise ValueError(f"need one goal box per environment ({self.n_envs}), got {ne}")
        rew = np.zeros(ne, np.float64)
        ins = np.zeros(ne, np.int64)
        call = lib().gg_goal_reward_noalloc if noalloc else lib().gg_goal_reward
        _check(call(self._h, bx.ctypes.data_as(C.c_void_p), rew.ctypes.data_as(C.c_void_p),
                    ins.ctypes.data_as(C.c_void_p), GG_MEM_HOST))
        return rew, ins

    def backward(self, dL_dx=None, dL_dv=None, n_steps=None):
        """Gradients of the last (differentiable) step call: returns
        (dL/dx0, dL/dv0, dL/dtwists) as NumPy arrays given dL/dx, dL/dv of the
        final state (None = zero)."""
        n = self.n
        gx = None if dL_dx is None else np.ascontiguousarray(dL_dx, np.float32).reshape(n, 3)
        gv = None if dL_dv is None else np.ascontiguousarray(dL_dv, np.float32).reshape(n, 3)
        ox = np.zeros((n, 3), np.float32)
        ov = np.zeros((n, 3), np.float32)
        steps = self.last_steps if n_steps is None else n_steps
        ot = np.zeros((steps, self.n_bodies, 6), np.float32)
        p = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
        _check(lib().gg_step_backward(self._h, p(gx), p(gv), p(ox), p(ov), p(ot) if ot.size else None,
                                      GG_MEM_HOST))
        return ox, ov, ot


def scene_sim(scene, **kw):
    """Sim initialised from a scenes.Scene (host arrays)."""
    args = dict(dt=scene.dt, alpha=scene.alpha, mu=scene.mu, n_iters=scene.n_iters,
                gravity=scene.gravity, env_offsets=scene.env_offsets)
    args.update(kw)
    return Sim(scene.x, scene.v, scene.radius, scene.bodies, **args)


def rollout_function():
    """torch.autograd.Function over a differentiable rollout:
    (x0, v0, twists) -> (x_final, v_final).  Each forward builds a simulation
    from (x0, v0) with GG_FLAG_TAPE, runs len(twists) steps and keeps it for the
    backward, which calls gg_step_backward (checkpointed recompute + adjoint
    kernels).  ``setup`` carries radius, bodies and Sim keyword arguments."""
    import torch

    class Rollout(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x0, v0, twists, setup):
            sim = Sim(x0.detach().cpu().numpy(), v0.detach().cpu().numpy(), setup["radius"], setup["bodies"],
                      differentiable=True, **setup.get("kwargs", {}))
            tw = twists.detach().cpu().numpy().astype(np.float32)
            sim.step(tw.shape[0], twists=tw)
            ctx.sim = sim
            x = torch.from_numpy(sim.read("pos")).to(x0.device)
            v = torch.from_numpy(sim.read("vel")).to(x0.device)
            return x, v

        @staticmethod
        def backward(ctx, gx, gv):
            sim = ctx.sim
            ox, ov, ot = sim.backward(None if gx is None else gx.detach().cpu().numpy(),
                                      None if gv is None else gv.detach().cpu().numpy())
            sim.close()
            dev = gx.device if gx is not None else gv.device
            return (torch.from_numpy(ox).to(dev), torch.from_numpy(ov).to(dev), torch.from_numpy(ot).to(dev), None)

    return Rollout
