"""Gym-style bulldozing environment around the simulator (arXiv 2306.01369,
Sec. III-A, "Bulldozing").

A batch of independent environments in one simulation (the batched form: one
particle segment and one set of bodies per environment).  Each environment is
a walled square arena holding a pile of grains, a goal box along the far side
and a bulldozer blade, a box body driven by a track steering model: the action
(a_lin, a_yaw) in [-1, 1]^2 sets the forward speed along the blade's heading
(v_max a_lin) and the yaw rate (yaw_max a_yaw) about the vertical through the
blade's centre.  One environment step runs `substeps` simulator steps of `dt`
(0.01 s by default, the coarse step the paper trains with), then observes each
environment through an ego camera (perspective, riding on the blade and
looking ahead of it) and a sky camera (orthographic, looking down on the whole
arena), both rendered on the device, plus the blade's planar pose (x, y, yaw);
the reward is the goal-box reward (100/n per grain inside the box, -d/n per
grain outside it at distance d).

The paper's arena, vehicle model, camera placement and control period are not
given; the values here are choices of this environment, stated in the
constructor's arguments.  The default pile is about four grains deep: at the
coarse 10 ms step, 20 projected-Jacobi sweeps cannot hold up much taller
stacks, which then sink into themselves (the collapse of tall stacks the paper
reports for this step size) until contacts exceed their capacity.  For the
same reason grains that the kinematic blade drives into the pile overlap
their neighbours deeply -- more neighbours than a sphere can touch without
overlap, and some sink into the floor -- so the contact capacity defaults to
64 per grain rather than the packing bound.
"""
from __future__ import annotations

import math

import numpy as np

from . import gg, scenes


class BulldozerEnv:
    """Batched bulldozing environment.

    reset() -> obs; step(actions (n_envs, 2)) -> (obs, reward (n_envs,),
    done (n_envs,), info).  obs = {"ego": (n_envs, H, W) depth, "sky":
    (n_envs, H, W) depth, "pose": (n_envs, 3) blade x, y (arena frame), yaw}.
    With device_obs=True the depth images are torch tensors on the device the
    simulation runs on (no host copy)."""

    def __init__(self, n_envs=4, n_particles=8192, seed=0, r=0.004, arena=0.7, pile=0.4, dt=0.01,
                 substeps=5, n_iters=20, mu=0.5, alpha=0.2, horizon=100, v_max=0.15, yaw_max=1.0,
                 blade=(0.015, 0.1, 0.05), ego=(64, 48), sky=(64, 64), ego_fov=70.0, graph=True,
                 precision=0, device_obs=False, max_contacts=64):
        self.n_envs, self.n_particles, self.r = int(n_envs), int(n_particles), float(r)
        self.arena, self.pile = float(arena), float(pile)
        self.dt, self.substeps, self.horizon = float(dt), int(substeps), int(horizon)
        self.v_max, self.yaw_max = float(v_max), float(yaw_max)
        self.blade = tuple(float(b) for b in blade)
        self.ego_size, self.sky_size, self.ego_fov = tuple(ego), tuple(sky), float(ego_fov)
        self.sim_kw = dict(dt=dt, n_iters=n_iters, mu=mu, alpha=alpha, graph=graph, precision=precision,
                           max_contacts=max_contacts)
        self.device_obs = bool(device_obs)
        self.seed = seed
        self.sim = None
        self._build(seed)

    # ---------------------------------------------------------------- layout
    def origin(self, e):
        """World position of environment e's arena corner (arenas on a grid,
        0.4 m apart)."""
        g = int(math.ceil(math.sqrt(self.n_envs)))
        pitch = self.arena + 0.4
        return (e % g) * pitch, (e // g) * pitch

    def goal_box(self, e):
        gx, gy = self.origin(e)
        a = self.arena
        return np.array([gx + 0.8 * a, gy, 0.0, gx + a, gy + a, 0.2], np.float32)

    def _build(self, seed):
        rng = np.random.default_rng(seed)
        xs, bodies, self.blade_index = [], [], []
        a, p = self.arena, self.pile
        for e in range(self.n_envs):
            gx, gy = self.origin(e)
            y0 = gy + 0.5 * (a - p)
            xs.append(scenes.packed_bed(self.n_particles, self.r, gx + 0.1 * a, gx + 0.1 * a + p, y0, y0 + p, rng))
            bodies += scenes.walled_box(gx, gx + a, gy, gy + a, env=e)
            self.blade_index.append(len(bodies))
            # the blade reaches 2 cm below the floor: no grain can be caught under
            # it, and a grain pressed into its face stays nearer that face than
            # the bottom face (whose normal would push it into the floor)
            bodies.append(scenes.box_tool((gx + 0.035, gy + 0.5 * a, self.blade[2] - 0.02), self.blade, env=e))
        self.x0 = np.ascontiguousarray(np.concatenate(xs), np.float32)
        self.radius = np.full(len(self.x0), self.r, np.float32)
        self.offsets = np.arange(self.n_envs + 1, dtype=np.int64) * self.n_particles
        self.bodies = bodies
        self.boxes = np.stack([self.goal_box(e) for e in range(self.n_envs)])
        # cameras: [ego_0, sky_0, ego_1, sky_1, ...]; the sky cameras never move
        cams = []
        for e in range(self.n_envs):
            gx, gy = self.origin(e)
            cams.append(scenes.perspective_camera((0, 0, 1), (1, 0, 1), self.ego_fov, self.ego_size[0],
                                                  self.ego_size[1], 1.0, env=e))
            cams.append(scenes.sky_camera(gx, gx + a, gy, gy + a, 0.4, self.sky_size[0], self.sky_size[1], env=e))
        self.cams = cams
        self.cam_array = gg.make_cameras(cams)
        self.cam_view = np.ctypeslib.as_array(self.cam_array)   # writes go to the camera array
        self.corners = np.array([self.origin(e) for e in range(self.n_envs)], np.float64)
        self.ego_px = self.ego_size[0] * self.ego_size[1]
        self.sky_px = self.sky_size[0] * self.sky_size[1]

    # ---------------------------------------------------------------- control
    def _ego_poses(self):
        """Ego camera poses (n_envs, 3, 4): 6 cm behind and 10 cm above the
        blade's top, looking at the floor 25 cm ahead of it."""
        x, y, th = self.state[:, 0], self.state[:, 1], self.state[:, 2]
        c, s = np.cos(th), np.sin(th)
        z = self.blade[2] - 0.02
        eye = np.stack([x - 0.06 * c, y - 0.06 * s, np.full_like(x, z + 0.10)], axis=1)
        tgt = np.stack([x + 0.25 * c, y + 0.25 * s, np.zeros_like(x)], axis=1)
        f = tgt - eye
        f /= np.linalg.norm(f, axis=1, keepdims=True)
        xa = np.cross(f, np.array([0.0, 0.0, 1.0]))
        xa /= np.linalg.norm(xa, axis=1, keepdims=True)
        ya = np.cross(f, xa)
        return np.concatenate([np.stack([xa, ya, f], axis=2), eye[:, :, None]], axis=2)

    def _twists(self, actions):
        """Per-substep body twists (substeps, n_bodies, 6) and the blade poses
        they lead to (the library advances t += dt nu, yaw += dt omega).  The
        vehicle stops where a step would bring the blade's centre closer to a
        wall than its half width plus 2 cm (it may still turn there, and move
        away from the wall), so the blade never crushes grains against the
        walls."""
        act = np.clip(np.asarray(actions, np.float64).reshape(self.n_envs, 2), -1.0, 1.0)
        tw = np.zeros((self.substeps, len(self.bodies), 6), np.float32)
        m = math.hypot(self.blade[0], self.blade[1]) + 0.02
        lo = self.corners + m
        hi = self.corners + self.arena - m

        def out(p):
            return (np.maximum(np.maximum(lo - p, p - hi), 0.0)).sum(axis=1)
        v0, w = self.v_max * act[:, 0], self.yaw_max * act[:, 1]
        b = np.asarray(self.blade_index)
        for k in range(self.substeps):
            xy, th = self.state[:, :2], self.state[:, 2]
            head = np.stack([np.cos(th), np.sin(th)], axis=1)
            v = np.where(out(xy + self.dt * v0[:, None] * head) > out(xy), 0.0, v0)
            nu = (v[:, None] * head).astype(np.float32)
            om = w.astype(np.float32)
            tw[k, b, 0:2] = nu
            tw[k, b, 5] = om
            self.state[:, 0:2] += self.dt * nu.astype(np.float64)
            self.state[:, 2] += self.dt * om.astype(np.float64)
        return tw

    # ---------------------------------------------------------------- Gym API
    def reset(self, seed=None):
        if seed is not None and seed != self.seed:
            self.seed = seed
            self._build(seed)
        if self.sim is not None:
            self.sim.close()
        self.sim = gg.Sim(self.x0, np.zeros_like(self.x0), self.radius, self.bodies, env_offsets=self.offsets,
                          **self.sim_kw)
        self.state = self.initial_state()
        self.t = 0
        return self.observe()

    def initial_state(self):
        """Blade (x, y, yaw) per environment at reset, x and y as the library
        holds them (binary32)."""
        t = np.array([self.bodies[b]["t"][:2] for b in self.blade_index], np.float32).astype(np.float64)
        return np.concatenate([t, np.zeros((self.n_envs, 1))], axis=1)

    def observe(self):
        self.cam_view["pose"][0::2] = self._ego_poses().reshape(self.n_envs, 12)
        total = self.n_envs * (self.ego_px + self.sky_px)
        per = self.ego_px + self.sky_px
        if self.device_obs:
            import torch
            buf = torch.empty(total, dtype=torch.float32, device="cuda")
            self.sim.render_cameras(self.cam_array, 2 * self.n_envs, buf)
            view = buf.view(self.n_envs, per)
        else:
            buf = np.empty(total, np.float32)
            self.sim.render_cameras(self.cam_array, 2 * self.n_envs, buf)
            view = buf.reshape(self.n_envs, per)
        ego = view[:, :self.ego_px].reshape(self.n_envs, self.ego_size[1], self.ego_size[0])
        sky = view[:, self.ego_px:].reshape(self.n_envs, self.sky_size[1], self.sky_size[0])
        # the blade's planar pose as the library advanced it
        P = self.sim.read("body_poses")[self.blade_index].astype(np.float64)
        pose = np.stack([P[:, 0, 3] - self.corners[:, 0], P[:, 1, 3] - self.corners[:, 1],
                         np.arctan2(P[:, 1, 0], P[:, 0, 0])], axis=1)
        return {"ego": ego, "sky": sky, "pose": pose}

    def step(self, actions):
        tw = self._twists(actions)
        self.sim.step(self.substeps, tw)
        self.t += 1
        obs = self.observe()
        reward, inside = self.sim.goal_reward(self.boxes)
        done = np.full(self.n_envs, self.t >= self.horizon)
        return obs, reward, done, {"inside": inside, "t": self.t}

    def cameras(self):
        """The camera dicts of the last observation (ego poses as rendered)."""
        out = []
        for k, c in enumerate(self.cams):
            A = self.cam_array[k]
            out.append(dict(c, pose=np.array(A.pose[:], np.float32).reshape(3, 4)))
        return out

    def close(self):
        if self.sim is not None:
            self.sim.close()
            self.sim = None
