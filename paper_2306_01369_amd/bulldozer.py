"""Gym-style bulldozing environment around the simulator (arXiv 2306.01369,
Sec. V-A, "Bulldozing").

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
constructor's arguments.
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

    def __init__(self, n_envs=4, n_particles=8192, seed=0, r=0.004, arena=0.6, pile=0.3, dt=0.01,
                 substeps=5, n_iters=20, mu=0.5, alpha=0.2, horizon=100, v_max=0.25, yaw_max=1.5,
                 blade=(0.015, 0.1, 0.04), ego=(64, 48), sky=(64, 64), ego_fov=70.0, graph=True,
                 precision=0, device_obs=False):
        self.n_envs, self.n_particles, self.r = int(n_envs), int(n_particles), float(r)
        self.arena, self.pile = float(arena), float(pile)
        self.dt, self.substeps, self.horizon = float(dt), int(substeps), int(horizon)
        self.v_max, self.yaw_max = float(v_max), float(yaw_max)
        self.blade = tuple(float(b) for b in blade)
        self.ego_size, self.sky_size, self.ego_fov = tuple(ego), tuple(sky), float(ego_fov)
        self.sim_kw = dict(dt=dt, n_iters=n_iters, mu=mu, alpha=alpha, graph=graph, precision=precision)
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
        return np.array([gx + 0.75 * a, gy, 0.0, gx + a, gy + a, 0.2], np.float32)

    def _build(self, seed):
        rng = np.random.default_rng(seed)
        xs, bodies, self.blade_index = [], [], []
        a, p = self.arena, self.pile
        for e in range(self.n_envs):
            gx, gy = self.origin(e)
            y0 = gy + 0.5 * (a - p)
            xs.append(scenes.packed_bed(self.n_particles, self.r, gx + 0.2 * a, gx + 0.2 * a + p, y0, y0 + p, rng))
            bodies += scenes.walled_box(gx, gx + a, gy, gy + a, env=e)
            self.blade_index.append(len(bodies))
            bodies.append(scenes.box_tool((gx + 0.06, gy + 0.5 * a, self.blade[2] + 0.002), self.blade, env=e))
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
        self.ego_px = self.ego_size[0] * self.ego_size[1]
        self.sky_px = self.sky_size[0] * self.sky_size[1]

    # ---------------------------------------------------------------- control
    def _ego_pose(self, e):
        x, y, th = self.state[e]
        c, s = math.cos(th), math.sin(th)
        z = self.blade[2] + 0.002
        eye = (x - 0.06 * c, y - 0.06 * s, z + 0.10)
        tgt = (x + 0.25 * c, y + 0.25 * s, 0.0)
        return scenes.camera_pose(eye, tgt)

    def _twists(self, actions):
        """Per-substep body twists (substeps, n_bodies, 6) and the blade poses
        they lead to (the library advances t += dt nu, yaw += dt omega)."""
        act = np.clip(np.asarray(actions, np.float64).reshape(self.n_envs, 2), -1.0, 1.0)
        tw = np.zeros((self.substeps, len(self.bodies), 6), np.float32)
        for k in range(self.substeps):
            for e in range(self.n_envs):
                x, y, th = self.state[e]
                v, w = self.v_max * act[e, 0], self.yaw_max * act[e, 1]
                nu = np.float32([v * math.cos(th), v * math.sin(th), 0.0])
                om = np.float32(w)
                b = self.blade_index[e]
                tw[k, b, 0:3] = nu
                tw[k, b, 5] = om
                self.state[e] = (x + self.dt * float(nu[0]), y + self.dt * float(nu[1]), th + self.dt * float(om))
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
        self.state = []
        for e in range(self.n_envs):
            t = self.bodies[self.blade_index[e]]["t"]
            self.state.append((float(np.float32(t[0])), float(np.float32(t[1])), 0.0))
        self.t = 0
        return self.observe()

    def observe(self):
        for e in range(self.n_envs):
            pose = np.asarray(self._ego_pose(e), np.float32).reshape(12)
            A = self.cam_array[2 * e]
            for q in range(12):
                A.pose[q] = float(pose[q])
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
        pose = np.array([(x - self.origin(e)[0], y - self.origin(e)[1], th)
                         for e, (x, y, th) in enumerate(self.state)])
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
