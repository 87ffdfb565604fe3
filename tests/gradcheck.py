"""Reference directional derivatives of a rollout (tests only).

The map (x0, v0, per-step twists) -> loss(x_N, v_N) is evaluated with the
FP64 oracle.  Two references: central differences along a direction with
every step's contact set held at that of the unperturbed run, and the
oracle's forward-mode (dual-number) step, exact along the direction with the
unperturbed run's decisions, the adjoint's own convention.  The differences
validate the dual numbers on smooth cases; at scale the dual numbers are the
reference, because central differences average across the non-smooth points
of the projection (unloaded contacts sit at the normal clamp)."""
import numpy as np

import oracle as O


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def box_sdf(p, center, half):
    q = np.abs(p - center) - half
    out = np.linalg.norm(np.maximum(q, 0.0), axis=1)
    ins = np.minimum(np.max(q, axis=1), 0.0)
    return out + ins


def box_sdf_grad(p, center, half):
    d = p - center
    s = np.where(d < 0, -1.0, 1.0)
    q = np.abs(d) - half
    m = np.maximum(q, 0.0)
    L = np.linalg.norm(m, axis=1)
    g = np.zeros_like(p)
    outside = L > 0
    g[outside] = s[outside] * m[outside] / L[outside, None]
    a = np.argmax(q, axis=1)
    ins = ~outside
    g[ins, a[ins]] = s[ins, a[ins]]
    return g


class TargetLoss:
    """L = sum_i sigmoid(-SDF_target(x_i)/width) + c . sum_i v_i"""

    def __init__(self, center, half, width=1e-3, vel_weight=(0.0, 0.0, 0.0)):
        self.center = np.asarray(center, float)
        self.half = np.asarray(half, float)
        self.width = width
        self.c = np.asarray(vel_weight, float)

    def __call__(self, x, v):
        return float(np.sum(sigmoid(-box_sdf(x, self.center, self.half) / self.width)) + np.sum(v @ self.c))

    def grads(self, x, v):
        z = -box_sdf(x, self.center, self.half) / self.width
        sg = sigmoid(z)
        dz = sg * (1 - sg) * (-1.0 / self.width)
        gx = dz[:, None] * box_sdf_grad(x, self.center, self.half)
        gv = np.broadcast_to(self.c, v.shape).copy()
        return gx, gv


def oracle_rollout(x0, v0, r, bodies, twists, detail=False, fixed=None, **kw):
    """Run the oracle; returns final state and, with detail, each step's
    (contact list, pair count).  fixed: such a list per step, held fixed."""
    orc = O.Oracle(x0, v0, r, bodies, **kw)
    lists = []
    for k in range(twists.shape[0]):
        orc.set_twists(twists[k], binary32=False)
        f = None if fixed is None else fixed[k]
        if detail or f is not None:
            d = orc.step(detail=True, fixed=f)
            lists.append((d["pairs"].copy(), d["n_pp"] if f is None else f[1]))
        else:
            orc.step()
    return orc.x, orc.v, lists


def fd_directional(loss, x0, v0, r, bodies, twists, d, h, **kw):
    """Central difference of loss along d with every step's contact set held at
    that of the unperturbed run (the adjoint's convention); also reports
    whether free detection would have kept the same sets."""
    dx, dv, dt = d
    x_, v_, base = oracle_rollout(x0, v0, r, bodies, twists, detail=True, **kw)
    xp, vp, _ = oracle_rollout(x0 + h * dx, v0 + h * dv, r, bodies, twists + h * dt, fixed=base, **kw)
    xm, vm, _ = oracle_rollout(x0 - h * dx, v0 - h * dv, r, bodies, twists - h * dt, fixed=base, **kw)
    _, _, free = oracle_rollout(x0 + h * dx, v0 + h * dv, r, bodies, twists + h * dt, detail=True, **kw)
    same = all(a[0].shape == b[0].shape and np.array_equal(a[0], b[0]) for a, b in zip(free, base))
    return (loss(xp, vp) - loss(xm, vm)) / (2 * h), same


def jvp_rollout(x0, v0, r, bodies, twists, dx0, dv0, dtwists, **kw):
    """Forward-mode rollout: final state and its tangent along (dx0, dv0,
    dtwists)."""
    orc = O.Oracle(x0, v0, r, bodies, **kw)
    orc.start_tangents(dx0, dv0)
    for k in range(twists.shape[0]):
        orc.set_twists(twists[k], binary32=False)
        orc.set_twist_tangents(dtwists[k])
        orc.step_jvp()
    return orc.x, orc.v, orc.dx, orc.dv


def jvp_directional(loss, x0, v0, r, bodies, twists, d, **kw):
    """Exact directional derivative of loss(x_N, v_N) along d = (dx, dv, dtw)."""
    dx, dv, dt = d
    xN, vN, dxN, dvN = jvp_rollout(x0, v0, r, bodies, twists, dx, dv, dt, **kw)
    gx, gv = loss.grads(xN, vN)
    return float(np.sum(gx * dxN) + np.sum(gv * dvN))
